"""Synthetic sparse-GLM instances with correlated Gaussian features.

Recipe (the paper's synthetic setting, Section 5.2; its generator sits in the
missing appendix, so the details below are this project's reading):

* rows of X are i.i.d. N(0, Sigma) with Sigma_ij = corr^|i-j|, drawn by the
  column recursion x_1 ~ N(0, 1), x_j = corr x_{j-1} + sqrt(1 - corr^2) e_j,
  which has exactly that covariance;
* each column is centred and scaled to unit population standard deviation
  (||x_j||^2 = n), then rounded to the storage type (f64, f32 or bf16 through
  f32), and every later quantity uses the rounded values;
* beta* has k_true entries equal to 1 at indices i * floor(p / k_true);
* noise is Gaussian with variance Var(X beta*) / SNR;
* least squares: y = X beta* + noise; logistic: y = sign(X beta* + noise) in
  {-1, +1} (sign 0 -> +1).

Draw order with ``numpy.random.default_rng(seed)``: all column innovations in
column order, then the noise.  X is stored column-major as a C-contiguous
``(p, n)`` array whose row j is column j.
"""
from dataclasses import dataclass, field
import math

import numpy as np


def round_bf16(a32: np.ndarray) -> np.ndarray:
    """float32 -> bf16 bit patterns (uint16), round to nearest even."""
    bits = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32)
    lsb = (bits >> np.uint32(16)) & np.uint32(1)
    r = (bits + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_to_f32(b16: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(b16, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


@dataclass
class Instance:
    name: str
    Xcm: np.ndarray          # (p, n) C-contiguous: column-major X in storage dtype
    y: np.ndarray            # (n,) float64
    n: int
    p: int
    loss: int                # 0 least squares, 1 logistic
    storage: str             # "f64" | "f32" | "bf16"
    beta_true: np.ndarray
    params: dict = field(default_factory=dict)

    def X64(self) -> np.ndarray:
        """Stored X exactly upcast to float64, column-major (p, n)."""
        if self.storage == "bf16":
            return bf16_to_f32(self.Xcm).astype(np.float64)
        return self.Xcm.astype(np.float64)


def make_instance(n, p, corr, k_true, snr, loss, seed, storage="f32", name="custom", **params):
    rng = np.random.default_rng(seed)
    if storage == "f64":
        Xcm = np.empty((p, n), dtype=np.float64)
    elif storage == "f32":
        Xcm = np.empty((p, n), dtype=np.float32)
    elif storage == "bf16":
        Xcm = np.empty((p, n), dtype=np.uint16)
    else:
        raise ValueError(storage)
    s = math.sqrt(1.0 - corr * corr)
    col = None
    for j in range(p):
        e = rng.standard_normal(n)
        col = e if col is None else corr * col + s * e
        c = col - col.mean()
        sd = c.std()
        c = c / sd if sd > 0 else c
        if storage == "f64":
            Xcm[j] = c
        elif storage == "f32":
            Xcm[j] = c.astype(np.float32)
        else:
            Xcm[j] = round_bf16(c.astype(np.float32))
    beta = np.zeros(p)
    step = p // k_true
    supp = [i * step for i in range(k_true)]
    beta[supp] = 1.0
    if storage == "bf16":
        cols = bf16_to_f32(Xcm[supp]).astype(np.float64)
    else:
        cols = Xcm[supp].astype(np.float64)
    signal = cols.sum(axis=0)
    sigma2 = signal.var() / snr
    noise = rng.standard_normal(n) * math.sqrt(sigma2)
    if loss == 0:
        y = signal + noise
    else:
        y = np.where(signal + noise >= 0.0, 1.0, -1.0)
    return Instance(name=name, Xcm=Xcm, y=np.ascontiguousarray(y, dtype=np.float64), n=n, p=p,
                    loss=loss, storage=storage, beta_true=beta, params=dict(params))


def make_nodes(p, m, seed, max_j0=64, max_j1=19):
    """m branch-and-bound nodes: |J0| ~ U{0..max_j0}, |J1| ~ U{0..max_j1},
    disjoint index sets drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    nodes = []
    for _ in range(m):
        n0 = int(rng.integers(0, max_j0 + 1))
        n1 = int(rng.integers(0, max_j1 + 1))
        idx = rng.choice(p, size=n0 + n1, replace=False)
        nodes.append((np.sort(idx[:n0]).astype(np.int32), np.sort(idx[n0:]).astype(np.int32)))
    return nodes


# Workloads: sizes, correlation, sparsity and loss of the measured configurations.
# M (box) is not stated for them; M = 2 is the paper's synthetic setting.
CONFIGS = {
    "ls_root_n500_p200_f64": dict(n=500, p=200, corr=0.5, k_true=10, snr=5.0, loss=0, seed=0,
                                  storage="f64", lambda2=1.0, k=10, M=2.0, tol=1e-8),
    "ls_root_n16384_p8192_f32": dict(n=16384, p=8192, corr=0.9, k_true=20, snr=5.0, loss=0, seed=0,
                                     storage="f32", lambda2=0.1, k=20, M=2.0, tol=1e-6),
    "logistic_root_n32768_p16384_f32": dict(n=32768, p=16384, corr=0.7, k_true=15, snr=5.0, loss=1,
                                            seed=0, storage="f32", lambda2=0.1, k=15, M=2.0,
                                            tol=1e-6),
    "ls_batch256_n16384_p8192_bf16": dict(n=16384, p=8192, corr=0.9, k_true=20, snr=5.0, loss=0,
                                          seed=0, storage="bf16", lambda2=0.1, k=20, M=2.0,
                                          tol=1e-6, m=256, node_seed=1),
}


def config_instance(name, **overrides):
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    keys = ("n", "p", "corr", "k_true", "snr", "loss", "seed", "storage")
    inst = make_instance(**{k: cfg[k] for k in keys}, name=name,
                         **{k: v for k, v in cfg.items() if k not in keys})
    return inst
