"""FP64 CPU oracle for the perspective-relaxation hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library never calls it, shares no code with it, and has no fallback to it.

All arrays are numpy float64 (vectors) plus the stored design matrix in its
storage dtype (column-major, i.e. a C-contiguous ``(p, n)`` array whose row j
is column j of X).  Function names follow the paper: ``g`` is g_N by Theorem compute_g_value,
``prox_gstar`` Algorithm 2, ``prox_g`` the Moreau identity (prox:gN), ``gstar``
the closed form of the conjugate, ``dual`` the Fenchel dual objective.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

FREE, ZERO, ONE = 0, 1, 2
LSQ, LOGISTIC = 0, 1
F64, F32, BF16 = 0, 1, 2
CONVERGED, MAXITER, INFEASIBLE, CUTOFF_PRUNE, CUTOFF_BRANCH = 1, 2, 3, 4, 5

_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_p = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_huber.restype = _d
        L.orc_huber.argtypes = [_d, _d]
        L.orc_prox_huber.restype = _d
        L.orc_prox_huber.argtypes = [_d, _d, _d]
        L.orc_g.restype = _d
        L.orc_g.argtypes = [_p, _p, _i64, _i32]
        L.orc_in_dom.restype = ctypes.c_int
        L.orc_in_dom.argtypes = [_p, _p, _i64, _i32, _d, _d]
        L.orc_gstar.restype = _d
        L.orc_gstar.argtypes = [_p, _p, _i64, _i32, _d]
        L.orc_prox_gstar.restype = None
        L.orc_prox_gstar.argtypes = [_p, _p, _i64, _d, _i32, _d, _p]
        L.orc_prox_g.restype = None
        L.orc_prox_g.argtypes = [_p, _p, _i64, _d, _i32, _d, _p]
        L.orc_loss.restype = _d
        L.orc_loss.argtypes = [ctypes.c_int, _p, _p, _i64]
        L.orc_loss_grad.restype = None
        L.orc_loss_grad.argtypes = [ctypes.c_int, _p, _p, _i64, _p]
        L.orc_neg_conj.restype = _d
        L.orc_neg_conj.argtypes = [ctypes.c_int, _p, _p, _i64]
        L.orc_matvec.restype = None
        L.orc_matvec.argtypes = [_p, ctypes.c_int, _i64, _i64, _p, _p]
        L.orc_rmatvec.restype = None
        L.orc_rmatvec.argtypes = [_p, ctypes.c_int, _i64, _i64, _p, _p]
        L.orc_power_norm2.restype = _d
        L.orc_power_norm2.argtypes = [_p, ctypes.c_int, _i64, _i64, _i64, _d]
        L.orc_primal.restype = _d
        L.orc_primal.argtypes = [_p, ctypes.c_int, _p, _i64, _i64, ctypes.c_int, _d, _d, _i32, _p, _p]
        L.orc_dual.restype = _d
        L.orc_dual.argtypes = [_p, ctypes.c_int, _p, _i64, _i64, ctypes.c_int, _d, _d, _i32, _p, _p]
        L.orc_solve.restype = ctypes.c_int
        L.orc_solve.argtypes = [_p, ctypes.c_int, _p, _i64, _i64, ctypes.c_int, _d, _d, _i32, _p,
                                _d, _d, _d, _i64, _d, _p, _p, _p, _p, _p, _i64, ctypes.c_int, _p, _p, _i64]
        L.orc_solve_acfgm.restype = ctypes.c_int
        L.orc_solve_acfgm.argtypes = [_p, ctypes.c_int, _p, _i64, _i64, ctypes.c_int, _d, _d, _i32, _p,
                                      _d, _d, _d, ctypes.c_int, _d, _d, _i64, _p, _p, _p, _p, _p, _p, _p, _p,
                                      _i64]
        L.orc_solve_bt.restype = ctypes.c_int
        L.orc_solve_bt.argtypes = [_p, ctypes.c_int, _p, _i64, _i64, ctypes.c_int, _d, _d, _i32, _p,
                                   _d, _d, _d, ctypes.c_int, _d, _d, _i64, _d, _p, _p, _p, _p, _p, _p, _p, _i64]
        L.orc_lasso_G.restype = _d
        L.orc_lasso_G.argtypes = [ctypes.c_int, _p, _i64, _d]
        L.orc_lasso_Gstar.restype = _d
        L.orc_lasso_Gstar.argtypes = [ctypes.c_int, _p, _i64, _d]
        L.orc_lasso_prox.restype = None
        L.orc_lasso_prox.argtypes = [ctypes.c_int, _p, _i64, _d, _d, _p]
        L.orc_lasso_dual.restype = _d
        L.orc_lasso_dual.argtypes = [_p, ctypes.c_int, _p, _i64, _i64, ctypes.c_int, _d, _p, _p]
        L.orc_lasso_solve.restype = ctypes.c_int
        L.orc_lasso_solve.argtypes = [_p, ctypes.c_int, _p, _i64, _i64, ctypes.c_int, _d, _d, _d, _d, _i64,
                                      ctypes.c_int, _p, _p, _p, _p, _p, _p, _i64]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _st(status, p):
    if status is None:
        return np.zeros(p, dtype=np.int8)
    s = np.ascontiguousarray(status, dtype=np.int8)
    assert s.shape == (p,)
    return s


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _xinfo(Xcm):
    """(pointer-holding array, dtype code, n, p) for a column-major matrix
    given as a C-contiguous (p, n) array (float64, float32 or uint16 bf16 bits)."""
    X = np.ascontiguousarray(Xcm)
    if X.dtype == np.float64:
        code = F64
    elif X.dtype == np.float32:
        code = F32
    elif X.dtype == np.uint16:
        code = BF16
    else:
        raise TypeError(f"unsupported matrix dtype {X.dtype}")
    p, n = X.shape
    return X, code, n, p


def status_vector(p, J0=(), J1=()):
    s = np.zeros(p, dtype=np.int8)
    s[list(J0)] = ZERO
    s[list(J1)] = ONE
    return s


def huber(a, M):
    return lib().orc_huber(float(a), float(M))


def prox_huber(u, c, M):
    return lib().orc_prox_huber(float(u), float(c), float(M))


def g(beta, k, status=None):
    b = _f64(beta)
    s = _st(status, b.size)
    return lib().orc_g(_ptr(b), _ptr(s), b.size, int(k))


def in_dom(beta, k, M, status=None, rtol=1e-9):
    b = _f64(beta)
    s = _st(status, b.size)
    return bool(lib().orc_in_dom(_ptr(b), _ptr(s), b.size, int(k), float(M), float(rtol)))


def gstar(alpha, k, M, status=None):
    a = _f64(alpha)
    s = _st(status, a.size)
    return lib().orc_gstar(_ptr(a), _ptr(s), a.size, int(k), float(M))


def prox_gstar(b, rho, k, M, status=None):
    b = _f64(b)
    s = _st(status, b.size)
    out = np.empty_like(b)
    lib().orc_prox_gstar(_ptr(b), _ptr(s), b.size, float(rho), int(k), float(M), _ptr(out))
    return out


def prox_g(v, rho, k, M, status=None):
    v = _f64(v)
    s = _st(status, v.size)
    out = np.empty_like(v)
    lib().orc_prox_g(_ptr(v), _ptr(s), v.size, float(rho), int(k), float(M), _ptr(out))
    return out


def loss(kind, u, y):
    u = _f64(u)
    y = _f64(y)
    return lib().orc_loss(int(kind), _ptr(u), _ptr(y), u.size)


def loss_grad(kind, u, y):
    u = _f64(u)
    y = _f64(y)
    out = np.empty_like(u)
    lib().orc_loss_grad(int(kind), _ptr(u), _ptr(y), u.size, _ptr(out))
    return out


def neg_conj(kind, zeta, y):
    z = _f64(zeta)
    y = _f64(y)
    return lib().orc_neg_conj(int(kind), _ptr(z), _ptr(y), z.size)


def matvec(Xcm, b):
    X, code, n, p = _xinfo(Xcm)
    b = _f64(b)
    out = np.empty(n)
    lib().orc_matvec(_ptr(X), code, n, p, _ptr(b), _ptr(out))
    return out


def rmatvec(Xcm, r):
    X, code, n, p = _xinfo(Xcm)
    r = _f64(r)
    out = np.empty(p)
    lib().orc_rmatvec(_ptr(X), code, n, p, _ptr(r), _ptr(out))
    return out


def power_norm2(Xcm, max_iter=2000, tol=1e-12):
    X, code, n, p = _xinfo(Xcm)
    return lib().orc_power_norm2(_ptr(X), code, n, p, int(max_iter), float(tol))


def primal(Xcm, y, beta, kind, lambda2, M, k, status=None):
    X, code, n, p = _xinfo(Xcm)
    y = _f64(y)
    b = _f64(beta)
    s = _st(status, p)
    return lib().orc_primal(_ptr(X), code, _ptr(y), n, p, int(kind), float(lambda2), float(M),
                            int(k), _ptr(s), _ptr(b))


def dual(Xcm, y, zeta, kind, lambda2, M, k, status=None):
    X, code, n, p = _xinfo(Xcm)
    y = _f64(y)
    z = _f64(zeta)
    s = _st(status, p)
    return lib().orc_dual(_ptr(X), code, _ptr(y), n, p, int(kind), float(lambda2), float(M),
                          int(k), _ptr(s), _ptr(z))


FISTA_GAP, FISTA, FISTA_FV, PGD = 0, 1, 2, 3


def solve(Xcm, y, kind, lambda2, M, k, status=None, L=0.0, tol=1e-8, eta=math.exp(3.0),
          max_iter=100000, cutoff=float("nan"), beta0=None, trace_cap=0, method=FISTA_GAP, restart_cap=0):
    """FISTA + duality-gap restart (or, with `method`, FISTA without restart,
    FISTA with function-value restart, or PGD).  Returns a dict with lb, ub,
    rel_gap, L, iters, restarts, status, beta, zeta (dual vector attaining
    lb), with trace_cap > 0 the traces of Phi - Psi and Phi per iterate, and
    with restart_cap > 0 the iterate indices at which restarts were taken."""
    X, code, n, p = _xinfo(Xcm)
    y = _f64(y)
    s = _st(status, p)
    b0 = None if beta0 is None else _f64(beta0)
    beta = np.empty(p)
    zeta = np.empty(n)
    res = np.zeros(8)
    trace = np.full(max(trace_cap, 1), np.nan)
    phi = np.full(max(trace_cap, 1), np.nan)
    rst = np.full(max(restart_cap, 1), -1, dtype=np.int64)
    lib().orc_solve(_ptr(X), code, _ptr(y), n, p, int(kind), float(lambda2), float(M), int(k),
                    _ptr(s), float(L), float(tol), float(eta), int(max_iter), float(cutoff),
                    None if b0 is None else _ptr(b0), _ptr(beta), _ptr(zeta), _ptr(res),
                    _ptr(trace) if trace_cap > 0 else None, int(trace_cap), int(method),
                    _ptr(phi) if trace_cap > 0 else None, _ptr(rst) if restart_cap > 0 else None,
                    int(restart_cap))
    m = int(res[4]) + 1
    return dict(lb=res[0], ub=res[1], rel_gap=res[2], L=res[3], iters=int(res[4]),
                restarts=int(res[5]), status=int(res[6]), beta=beta, zeta=zeta,
                trace=trace[:m] if trace_cap > 0 else None, phi_trace=phi[:m] if trace_cap > 0 else None,
                restart_at=rst[:min(int(res[5]), restart_cap)] if restart_cap > 0 else None)


def num_threads():
    return lib().orc_num_threads()


def solve_acfgm(Xcm, y, kind, lambda2, M, k, status=None, L0=1.0, c=2.0, b=0.1, restart=True, tol=1e-8,
                eta=math.exp(3.0), max_iter=100000, beta0=None, trace_cap=0):
    """AC-FGM (Li and Lan) with, if `restart`, the duality-gap restart.
    Returns lb, ub, rel_gap, L1 (accepted first-step constant), iters
    (evaluations), restarts, status, rejected (line-search trials), beta (the
    iterate attaining ub), zeta (dual vector attaining lb), and with
    trace_cap > 0 per-evaluation traces: gap, phi, lhat, step (epoch step
    index t, negative for a rejected trial)."""
    X, code, n, p = _xinfo(Xcm)
    y = _f64(y)
    s = _st(status, p)
    b0 = None if beta0 is None else _f64(beta0)
    beta = np.empty(p)
    zeta = np.empty(n)
    res = np.zeros(8)
    tr = [np.full(max(trace_cap, 1), np.nan) for _ in range(4)]
    lib().orc_solve_acfgm(_ptr(X), code, _ptr(y), n, p, int(kind), float(lambda2), float(M), int(k), _ptr(s),
                          float(L0), float(c), float(b), int(bool(restart)), float(tol), float(eta), int(max_iter),
                          None if b0 is None else _ptr(b0), _ptr(beta), _ptr(zeta), _ptr(res),
                          *[(_ptr(a) if trace_cap > 0 else None) for a in tr], int(trace_cap))
    m = int(res[4]) + 1
    out = dict(lb=res[0], ub=res[1], rel_gap=res[2], L1=res[3], iters=int(res[4]), restarts=int(res[5]),
               status=int(res[6]), rejected=int(res[7]), beta=beta, zeta=zeta)
    if trace_cap > 0:
        out.update(trace=tr[0][:m], phi_trace=tr[1][:m], lhat=tr[2][:m], step=tr[3][:m])
    return out


def solve_bt(Xcm, y, kind, lambda2, M, k, status=None, L0=1.0, c=2.0, Lmax=None, restart=True, tol=1e-8,
             eta=math.exp(3.0), max_iter=100000, cutoff=float("nan"), beta0=None, trace_cap=0):
    """FISTA with backtracking (Beck's monotone rule from L0, factor c, capped
    at Lmax: default the loss curvature times ||X||_2^2 by power iteration)
    and, if `restart`, the duality-gap restart.  Returns lb, ub, rel_gap, L
    (final), iters (accepted), restarts, status, rejected, beta (last
    iterate), zeta (dual vector attaining lb), and with trace_cap > 0 per
    accepted iterate: trace (gap), phi_trace, L_trace."""
    X, code, n, p = _xinfo(Xcm)
    y = _f64(y)
    s = _st(status, p)
    if Lmax is None:
        nrm = lib().orc_power_norm2(_ptr(X), code, n, p, 2000, 1e-12)
        Lmax = (2.0 if kind == LSQ else 0.25) * nrm
    b0 = None if beta0 is None else _f64(beta0)
    beta = np.empty(p)
    zeta = np.empty(n)
    res = np.zeros(8)
    tr = [np.full(max(trace_cap, 1), np.nan) for _ in range(3)]
    rc = lib().orc_solve_bt(_ptr(X), code, _ptr(y), n, p, int(kind), float(lambda2), float(M), int(k), _ptr(s),
                            float(L0), float(c), float(Lmax), int(bool(restart)), float(tol), float(eta),
                            int(max_iter), float(cutoff), None if b0 is None else _ptr(b0), _ptr(beta), _ptr(zeta),
                            _ptr(res), *[(_ptr(a) if trace_cap > 0 else None) for a in tr], int(trace_cap))
    if rc < 0:
        raise ValueError("solve_bt: needs L0 > 0, c > 1 and Lmax >= L0")
    m = int(res[4]) + 1
    out = dict(lb=res[0], ub=res[1], rel_gap=res[2], L=res[3], iters=int(res[4]), restarts=int(res[5]),
               status=int(res[6]), rejected=int(res[7]), beta=beta, zeta=zeta, Lmax=float(Lmax))
    if trace_cap > 0:
        out.update(trace=tr[0][:m], phi_trace=tr[1][:m], L_trace=tr[2][:m])
    return out


L1_REG, L1_BALL = 0, 1


def lasso_G(kind, beta, lam):
    b = _f64(beta)
    return lib().orc_lasso_G(int(kind), _ptr(b), b.size, float(lam))


def lasso_Gstar(kind, w, lam):
    a = _f64(w)
    return lib().orc_lasso_Gstar(int(kind), _ptr(a), a.size, float(lam))


def lasso_prox(kind, v, t, lam):
    v = _f64(v)
    out = np.empty_like(v)
    lib().orc_lasso_prox(int(kind), _ptr(v), v.size, float(t), float(lam), _ptr(out))
    return out


def lasso_dual(Xcm, y, kind, lam, zeta):
    """(Psi, scale) at the dual-feasible point built from zeta (see oracle.c)."""
    X, code, n, p = _xinfo(Xcm)
    y = _f64(y)
    z = _f64(zeta)
    sc = np.zeros(1)
    v = lib().orc_lasso_dual(_ptr(X), code, _ptr(y), n, p, int(kind), float(lam), _ptr(z), _ptr(sc))
    return v, float(sc[0])


def lasso_solve(Xcm, y, kind, lam, L=0.0, tol=1e-8, eta=math.exp(3.0), max_iter=100000, method=FISTA_GAP,
                beta0=None, trace_cap=0):
    """FISTA (with the duality-gap restart unless method == FISTA) on the LASSO
    problem of `kind` (L1_REG: ||y - X b||^2 + lam ||b||_1; L1_BALL: the same
    loss over ||b||_1 <= lam).  Returns lb, ub, rel_gap, L, iters, restarts,
    status, beta (iterate attaining ub), zeta (dual point attaining lb),
    traces of gap and Phi with trace_cap > 0."""
    X, code, n, p = _xinfo(Xcm)
    y = _f64(y)
    b0 = None if beta0 is None else _f64(beta0)
    beta = np.empty(p)
    zeta = np.empty(n)
    res = np.zeros(8)
    trace = np.full(max(trace_cap, 1), np.nan)
    phi = np.full(max(trace_cap, 1), np.nan)
    lib().orc_lasso_solve(_ptr(X), code, _ptr(y), n, p, int(kind), float(lam), float(L), float(tol), float(eta),
                          int(max_iter), int(method), None if b0 is None else _ptr(b0), _ptr(beta), _ptr(zeta),
                          _ptr(res), _ptr(trace) if trace_cap > 0 else None,
                          _ptr(phi) if trace_cap > 0 else None, int(trace_cap))
    m = int(res[4]) + 1
    return dict(lb=res[0], ub=res[1], rel_gap=res[2], L=res[3], iters=int(res[4]), restarts=int(res[5]),
                status=int(res[6]), beta=beta, zeta=zeta,
                trace=trace[:m] if trace_cap > 0 else None, phi_trace=phi[:m] if trace_cap > 0 else None)
