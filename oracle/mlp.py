"""FP64 CPU oracle for the learned warm start (per-coordinate MLP).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may use it; the product library shares
no code with it and never calls it.

The learned part is not in the paper: it proposes a starting point for a
child node of branch and bound from its parent's solution, and the solver's
FP64 duality gap decides whether that start is used, so no bound depends on
it.  Everything here is plain numpy in float64, written from the definitions:

* features of coordinate j of a child node, from the parent solution beta and
  h = X^T (y - X beta) (least squares):
      f0 = beta_j
      f1 = h_j / max_i |h_i|            (0 if h = 0)
      f2 = #{i : |beta_i| > |beta_j|} / p
      f3 = child status of j: -1 fixed to zero, 0 free, +1 fixed to one
      f4 = lambda2
      f5 = |J1| / k,  f6 = |J0| / k,  f7 = kbar / k,  kbar = min(k - |J1|, #free)
* network 8 -> 64 -> 64 -> 1 with ReLU, flat parameter vector
      W1 (64 x 8) | b1 (64) | W2 (64 x 64) | b2 (64) | w3 (64) | b3 (1)   = 4801
  (row-major weights, out = w3 . relu(W2 relu(W1 f + b1) + b2) + b3);
* the network predicts the change of each coordinate from parent to child;
  loss = mean over rows of (out - t)^2, t = beta_child_j - beta_parent_j;
* Adam (Kingma and Ba 2015) with bias correction.
"""
import numpy as np

NF, H = 8, 64
OFF_W1, OFF_B1 = 0, 512
OFF_W2, OFF_B2 = 576, 4672
OFF_W3, OFF_B3 = 4736, 4800
NPARAM = 4801


def unpack(params):
    """Views (W1, b1, W2, b2, w3, b3) of a flat parameter vector."""
    P = np.asarray(params, dtype=np.float64)
    assert P.shape == (NPARAM,)
    return (P[OFF_W1:OFF_B1].reshape(H, NF), P[OFF_B1:OFF_W2], P[OFF_W2:OFF_B2].reshape(H, H),
            P[OFF_B2:OFF_W3], P[OFF_W3:OFF_B3], P[OFF_B3])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def forward(params, F):
    """Network output for every row of F (rows x 8)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    F = np.asarray(F, dtype=np.float64)
    a1 = np.maximum(F @ W1.T + b1, 0.0)
    a2 = np.maximum(a1 @ W2.T + b2, 0.0)
    return a2 @ w3 + b3


def loss_grad(params, F, T):
    """(loss, gradient) of loss = mean_r (out_r - T_r)^2 by backpropagation,
    each step the chain rule applied to one layer of forward()."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    F = np.asarray(F, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    N = F.shape[0]
    z1 = F @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    out = a2 @ w3 + b3
    d = out - T
    loss = float(np.mean(d * d)) if N else 0.0
    dout = 2.0 * d / max(N, 1)               # d loss / d out
    g_w3 = a2.T @ dout
    g_b3 = dout.sum()
    dz2 = np.outer(dout, w3) * (z2 > 0)      # d loss / d z2
    g_W2 = dz2.T @ a1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g_W1 = dz1.T @ F
    g_b1 = dz1.sum(axis=0)
    return loss, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (params, m, v)."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def features(beta, h, status, lambda2, k):
    """Feature rows (p x 8) of a child node; status uses the oracle's codes
    (0 free, 1 fixed to zero, 2 fixed to one)."""
    beta = np.asarray(beta, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    st = np.asarray(status)
    p = beta.size
    n0 = int(np.sum(st == 1))
    n1 = int(np.sum(st == 2))
    kbar = min(k - n1, int(np.sum(st == 0)))
    a = np.abs(beta)
    hmax = np.max(np.abs(h)) if p else 0.0
    F = np.zeros((p, NF))
    F[:, 0] = beta
    F[:, 1] = h / hmax if hmax > 0 else 0.0
    srt = np.sort(a)
    F[:, 2] = (p - np.searchsorted(srt, a, side="right")) / p   # count of strictly larger
    F[:, 3] = np.where(st == 1, -1.0, np.where(st == 2, 1.0, 0.0))
    F[:, 4] = lambda2
    F[:, 5] = n1 / k
    F[:, 6] = n0 / k
    F[:, 7] = kbar / k
    return F


def init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, NF)) * np.sqrt(6.0 / NF)
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    w3 = rng.uniform(-1, 1, H) * np.sqrt(6.0 / H) * 0.1
    return pack(W1, np.zeros(H), W2, np.zeros(H), w3, 0.0)
