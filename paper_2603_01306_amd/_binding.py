"""ctypes binding of libpr (include/pr.h).  Argument marshalling only: every
step of the solve runs in the HIP kernels of libpr.so.  torch is used for
device memory and the current stream.  Importing this module does not need a
GPU; calling into the library does, and there is no fallback when libpr.so
is missing."""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpr.so")

PR_OK, PR_EINVAL, PR_EOVERLAP, PR_EDEVICE, PR_ENOMEM = 0, -1, -2, -3, -4
PROX_NOALLOC_MAX_P = 1048576
DEBUG_GRAM_RECHECK, DEBUG_FORCE_BATCH = 1, 2
CONVERGED, MAXITER, INFEASIBLE, CUTOFF_PRUNE, CUTOFF_BRANCH = 1, 2, 3, 4, 5
FREE, ZERO, ONE = 0, 1, 2
FISTA_GAP, FISTA, FISTA_FV, PGD, ACFGM_GAP, ACFGM, FISTA_BT_GAP, FISTA_BT = 0, 1, 2, 3, 4, 5, 6, 7
L1_REG, L1_BALL = 0, 1
BNB_OPTIMAL, BNB_NODE_LIMIT, BNB_TIME_LIMIT = 1, 2, 3
LSQ, LOGISTIC = 0, 1
F64, F32, BF16 = 0, 1, 2

EXPORTS = ["pr_opts_default", "pr_ctx_create", "pr_ctx_destroy", "pr_ctx_norm2", "pr_ctx_enable_gram", "pr_solve",
           "pr_prox", "pr_regularizer", "pr_dual_bound", "pr_gemv", "pr_gemv_t", "pr_gemv_t2", "pr_solve_batch",
           "pr_time_gemv_t", "pr_time_gemv", "pr_time_read", "pr_time_batch_gemm", "pr_time_gram_gemm", "pr_batch_union_size", "pr_time_prox", "pr_batch_tuning", "pr_gemm", "pr_mlp_features", "pr_mlp_forward",
           "pr_mlp_workspace", "pr_mlp_grad", "pr_mlp_adam", "pr_mlp_warm_start", "pr_bnb_opts_default", "pr_bnb", "pr_prox_noalloc", "pr_ctx_set_debug", "pr_lasso_solve", "pr_strerror"]

MLP_NFEAT, MLP_NPARAM = 8, 4801


class PrProblem(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("xdtype", ctypes.c_int32), ("loss", ctypes.c_int32),
                ("y", ctypes.c_void_p), ("n", ctypes.c_int64), ("p", ctypes.c_int64)]


class PrNode(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("pad0", ctypes.c_int32), ("lambda2", ctypes.c_double),
                ("M", ctypes.c_double), ("J0", ctypes.c_void_p), ("n0", ctypes.c_int64),
                ("J1", ctypes.c_void_p), ("n1", ctypes.c_int64)]


class PrOpts(ctypes.Structure):
    _fields_ = [("rel_gap_tol", ctypes.c_double), ("eta", ctypes.c_double),
                ("cutoff", ctypes.c_double), ("L", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("method", ctypes.c_int32), ("pad0", ctypes.c_int32), ("trace", ctypes.c_void_p),
                ("acfgm_b", ctypes.c_double), ("acfgm_c", ctypes.c_double), ("L0", ctypes.c_double)]


class PrLasso(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad0", ctypes.c_int32), ("lam", ctypes.c_double)]


class PrBnbOpts(ctypes.Structure):
    _fields_ = [("rel_gap_tol", ctypes.c_double), ("time_limit_s", ctypes.c_double), ("max_nodes", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("node_opts", PrOpts)]


class PrBnbResult(ctypes.Structure):
    _fields_ = [("lower_bound", ctypes.c_double), ("upper_bound", ctypes.c_double), ("rel_gap", ctypes.c_double),
                ("seconds", ctypes.c_double), ("relaxation_seconds", ctypes.c_double),
                ("nodes_solved", ctypes.c_int64), ("nodes_pruned", ctypes.c_int64), ("nodes_open", ctypes.c_int64),
                ("max_depth", ctypes.c_int32), ("status", ctypes.c_int32)]


class PrResult(ctypes.Structure):
    _fields_ = [("lower_bound", ctypes.c_double), ("primal", ctypes.c_double),
                ("rel_gap", ctypes.c_double), ("L", ctypes.c_double), ("iters", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("status", ctypes.c_int32), ("trials", ctypes.c_int32)]

    def as_dict(self):
        return dict(lower_bound=self.lower_bound, primal=self.primal, rel_gap=self.rel_gap, L=self.L,
                    iters=self.iters, restarts=self.restarts, status=self.status, trials=self.trials)


_lib = None


def load():
    """Load libpr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libpr.so not found at {LIB_PATH}: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.pr_opts_default.restype = None
        L.pr_opts_default.argtypes = [ctypes.POINTER(PrOpts)]
        L.pr_ctx_create.restype = ctypes.c_int
        L.pr_ctx_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(PrProblem), ctypes.c_int32, P]
        L.pr_ctx_destroy.restype = ctypes.c_int
        L.pr_ctx_destroy.argtypes = [P]
        L.pr_ctx_set_debug.restype = ctypes.c_int
        L.pr_ctx_set_debug.argtypes = [P, ctypes.c_int32]
        L.pr_ctx_norm2.restype = ctypes.c_int
        L.pr_ctx_norm2.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
        L.pr_solve.restype = ctypes.c_int
        L.pr_solve.argtypes = [P, ctypes.POINTER(PrNode), ctypes.POINTER(PrOpts), P, P, P,
                               ctypes.POINTER(PrResult)]
        L.pr_prox.restype = ctypes.c_int
        L.pr_prox.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                              P, P]
        L.pr_prox_noalloc.restype = ctypes.c_int
        L.pr_prox_noalloc.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                      P, P]
        L.pr_regularizer.restype = ctypes.c_int
        L.pr_regularizer.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.pr_dual_bound.restype = ctypes.c_int
        L.pr_dual_bound.argtypes = [P, ctypes.POINTER(PrNode), P, P, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        L.pr_gemv.restype = ctypes.c_int
        L.pr_gemv.argtypes = [P, P, P]
        L.pr_gemv_t.restype = ctypes.c_int
        L.pr_gemv_t.argtypes = [P, P, P]
        L.pr_gemv_t2.restype = ctypes.c_int
        L.pr_gemv_t2.argtypes = [P, P, P, P, P]
        L.pr_time_gemv_t.restype = ctypes.c_int
        L.pr_time_gemv_t.argtypes = [P, P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.pr_time_gemv.restype = ctypes.c_int
        L.pr_time_gemv.argtypes = [P, P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.pr_time_read.restype = ctypes.c_int
        L.pr_time_read.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P,
                                   ctypes.POINTER(ctypes.c_double)]
        L.pr_lasso_solve.restype = ctypes.c_int
        L.pr_lasso_solve.argtypes = [P, ctypes.POINTER(PrLasso), ctypes.POINTER(PrOpts), P, P, P,
                                     ctypes.POINTER(PrResult)]
        L.pr_solve_batch.restype = ctypes.c_int
        L.pr_solve_batch.argtypes = [P, ctypes.POINTER(PrNode), ctypes.c_int32, ctypes.POINTER(PrOpts),
                                     P, P, ctypes.POINTER(PrResult)]
        L.pr_time_prox.restype = ctypes.c_int
        L.pr_time_prox.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double, P, P,
                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.pr_batch_tuning.restype = ctypes.c_int
        L.pr_batch_tuning.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.pr_time_batch_gemm.restype = ctypes.c_int
        L.pr_time_batch_gemm.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        L.pr_time_gram_gemm.restype = ctypes.c_int
        L.pr_time_gram_gemm.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.pr_batch_union_size.restype = ctypes.c_int
        L.pr_batch_union_size.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]
        L.pr_gemm.restype = ctypes.c_int
        L.pr_gemm.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_int32]
        L.pr_mlp_features.restype = ctypes.c_int
        L.pr_mlp_features.argtypes = [P, ctypes.POINTER(PrNode), ctypes.c_int32, P, P, P, P]
        L.pr_mlp_forward.restype = ctypes.c_int
        L.pr_mlp_forward.argtypes = [P, P, P, ctypes.c_int64, P]
        L.pr_mlp_workspace.restype = ctypes.c_int64
        L.pr_mlp_workspace.argtypes = [ctypes.c_int64]
        L.pr_mlp_grad.restype = ctypes.c_int
        L.pr_mlp_grad.argtypes = [P, P, P, P, ctypes.c_int64, P, P]
        L.pr_mlp_adam.restype = ctypes.c_int
        L.pr_mlp_adam.argtypes = [P, P, P, P, P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double]
        L.pr_mlp_warm_start.restype = ctypes.c_int
        L.pr_mlp_warm_start.argtypes = [P, ctypes.POINTER(PrNode), ctypes.c_int32, P, P, P,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
        L.pr_ctx_enable_gram.restype = ctypes.c_int
        L.pr_ctx_enable_gram.argtypes = [P]
        L.pr_bnb_opts_default.restype = None
        L.pr_bnb_opts_default.argtypes = [ctypes.POINTER(PrBnbOpts)]
        L.pr_bnb.restype = ctypes.c_int
        L.pr_bnb.argtypes = [P, ctypes.POINTER(PrNode), ctypes.POINTER(PrBnbOpts), P, ctypes.POINTER(PrBnbResult)]
        L.pr_strerror.restype = ctypes.c_char_p
        L.pr_strerror.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


class PrError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {load().pr_strerror(code).decode()} ({code})")
        self.code = code


def _check(code, what):
    if code != PR_OK:
        raise PrError(code, what)


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def default_opts(**kw):
    o = PrOpts()
    load().pr_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if v is None:
            continue
        if k == "trace":
            v = v.data_ptr()  # a float64 CUDA tensor of 2 * (max_iter + 1) entries
        setattr(o, k, v)
    return o


class Node:
    """A branch-and-bound node (k, lambda2, M, J0, J1); index arrays are kept alive here."""

    def __init__(self, k, lambda2, M=2.0, J0=(), J1=()):
        self.k = int(k)
        self.lambda2 = float(lambda2)
        self.M = float(M)
        self.J0 = np.ascontiguousarray(np.asarray(J0, dtype=np.int32).ravel())
        self.J1 = np.ascontiguousarray(np.asarray(J1, dtype=np.int32).ravel())

    def c(self):
        s = PrNode()
        s.k = self.k
        s.lambda2 = self.lambda2
        s.M = self.M
        s.J0 = self.J0.ctypes.data if self.J0.size else None
        s.n0 = self.J0.size
        s.J1 = self.J1.ctypes.data if self.J1.size else None
        s.n1 = self.J1.size
        return s

    def status(self, p):
        st = np.zeros(p, dtype=np.int8)
        st[self.J0] = ZERO
        st[self.J1] = ONE
        return st


def _xdtype(X):
    import torch
    if X.dtype == torch.float64:
        return F64
    if X.dtype == torch.float32:
        return F32
    if X.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported X dtype {X.dtype}")


class Context:
    """pr_ctx over a device-resident problem.  Xcm: CUDA tensor of shape (p, n)
    (row j = column j of X, i.e. column-major X), float64 / float32 / bfloat16;
    y: CUDA float64 tensor (n,)."""

    def __init__(self, Xcm, y, loss, max_batch=1):
        import torch
        assert Xcm.is_cuda and y.is_cuda and Xcm.is_contiguous() and y.is_contiguous()
        assert y.dtype == torch.float64
        self.X = Xcm
        self.y = y
        self.p, self.n = Xcm.shape
        self.loss = int(loss)
        self.max_batch = int(max_batch)
        prob = PrProblem()
        prob.X = Xcm.data_ptr()
        prob.xdtype = _xdtype(Xcm)
        prob.loss = self.loss
        prob.y = y.data_ptr()
        prob.n = self.n
        prob.p = self.p
        h = ctypes.c_void_p()
        _check(load().pr_ctx_create(ctypes.byref(h), ctypes.byref(prob), int(max_batch), _stream_ptr()),
               "pr_ctx_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().pr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def enable_gram(self):
        """Switch the context's least-squares solves to the Gram form h = b - G x."""
        _check(load().pr_ctx_enable_gram(self.h), "pr_ctx_enable_gram")

    def set_debug(self, flags):
        """Test switches (pr_ctx_set_debug); DEBUG_GRAM_RECHECK forces Gram-mode
        solves onto the matrix-vector re-solve."""
        _check(load().pr_ctx_set_debug(self.h, int(flags)), "pr_ctx_set_debug")

    def norm2(self):
        v = ctypes.c_double()
        _check(load().pr_ctx_norm2(self.h, ctypes.byref(v)), "pr_ctx_norm2")
        return v.value

    def solve(self, node, beta0=None, want_beta=True, want_zeta=False, **opts):
        import torch
        o = default_opts(**opts)
        dev = self.X.device
        beta = torch.empty(self.p, dtype=torch.float64, device=dev) if want_beta else None
        zeta = torch.empty(self.n, dtype=torch.float64, device=dev) if want_zeta else None
        if beta0 is not None:
            beta0 = beta0.to(device=dev, dtype=torch.float64).contiguous()
        res = PrResult()
        nd = node.c()
        _check(load().pr_solve(self.h, ctypes.byref(nd), ctypes.byref(o), _dptr(beta0), _dptr(beta),
                               _dptr(zeta), ctypes.byref(res)), "pr_solve")
        out = res.as_dict()
        out["beta"] = beta
        out["zeta"] = zeta
        return out

    def lasso_solve(self, kind, lam, beta0=None, want_beta=True, want_zeta=False, **opts):
        """LASSO with the duality-gap restart (kind L1_REG: penalty lam; L1_BALL:
        radius lam) on the context's least-squares problem."""
        import torch
        o = default_opts(**opts)
        dev = self.X.device
        beta = torch.empty(self.p, dtype=torch.float64, device=dev) if want_beta else None
        zeta = torch.empty(self.n, dtype=torch.float64, device=dev) if want_zeta else None
        if beta0 is not None:
            beta0 = beta0.to(device=dev, dtype=torch.float64).contiguous()
        lp = PrLasso()
        lp.kind = int(kind)
        lp.lam = float(lam)
        res = PrResult()
        _check(load().pr_lasso_solve(self.h, ctypes.byref(lp), ctypes.byref(o), _dptr(beta0), _dptr(beta),
                                     _dptr(zeta), ctypes.byref(res)), "pr_lasso_solve")
        out = res.as_dict()
        out["beta"] = beta
        out["zeta"] = zeta
        return out

    def solve_batch(self, nodes, B0=None, want_beta=True, **opts):
        import torch
        o = default_opts(**opts)
        m = len(nodes)
        arr = (PrNode * m)(*[nd.c() for nd in nodes])
        res = (PrResult * m)()
        dev = self.X.device
        Bout = torch.empty((m, self.p), dtype=torch.float64, device=dev) if want_beta else None
        if B0 is not None:
            B0 = B0.to(device=dev, dtype=torch.float64).contiguous()
        _check(load().pr_solve_batch(self.h, arr, m, ctypes.byref(o), _dptr(B0), _dptr(Bout), res),
               "pr_solve_batch")
        return [r.as_dict() for r in res], Bout

    def batch_tuning(self, tiles):
        """Autotuned (forward, transpose) split counts for 1 .. tiles active 64-row tiles."""
        a = (ctypes.c_int32 * tiles)()
        b = (ctypes.c_int32 * tiles)()
        _check(load().pr_batch_tuning(self.h, int(tiles), a, b), "pr_batch_tuning")
        return list(a), list(b)

    def time_batch_gemm(self, m, reps=20):
        """(ms forward GEMM, ms transpose GEMM) per launch for a batch of m nodes."""
        a = ctypes.c_double()
        b = ctypes.c_double()
        _check(load().pr_time_batch_gemm(self.h, int(m), int(reps), ctypes.byref(a), ctypes.byref(b)),
               "pr_time_batch_gemm")
        return a.value, b.value

    def time_gram_gemm(self, m, reps=20):
        """ms per launch of the batched Gram product G X_it for m active nodes."""
        a = ctypes.c_double()
        _check(load().pr_time_gram_gemm(self.h, int(m), int(reps), ctypes.byref(a)), "pr_time_gram_gemm")
        return a.value

    def batch_union_size(self):
        """(|U|, padded size, nonzeros outside U at the nodes' last iterates)
        of the support union the last batched Gram solve compacted its product
        to, (0, 0, 0) when it ran without."""
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        o = ctypes.c_int64()
        _check(load().pr_batch_union_size(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(o)),
               "pr_batch_union_size")
        return a.value, b.value, o.value

    def bnb(self, root, node_opts=None, **opts):
        """Branch and bound from `root`; returns (result dict, incumbent (p,) float64)."""
        import torch
        o = PrBnbOpts()
        load().pr_bnb_opts_default(ctypes.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        if node_opts:
            o.node_opts = default_opts(**node_opts)
        beta = torch.zeros(self.p, dtype=torch.float64, device=self.X.device)
        res = PrBnbResult()
        nd = root.c()
        _check(load().pr_bnb(self.h, ctypes.byref(nd), ctypes.byref(o), _dptr(beta), ctypes.byref(res)), "pr_bnb")
        out = {f: getattr(res, f) for f, _ in PrBnbResult._fields_}
        return out, beta

    def mlp_features(self, nodes, Bparent, Bchild=None):
        """Feature rows (m*p, 8) bfloat16 of child nodes from their parents'
        solutions (m, p) float64; with Bchild also the targets (m*p,) float32."""
        import torch
        m = len(nodes)
        dev = self.X.device
        arr = (PrNode * m)(*[nd.c() for nd in nodes])
        Bparent = Bparent.to(device=dev, dtype=torch.float64).contiguous()
        F = torch.empty((m * self.p, MLP_NFEAT), dtype=torch.bfloat16, device=dev)
        T = None
        if Bchild is not None:
            Bchild = Bchild.to(device=dev, dtype=torch.float64).contiguous()
            T = torch.empty(m * self.p, dtype=torch.float32, device=dev)
        _check(load().pr_mlp_features(self.h, arr, m, _dptr(Bparent), _dptr(Bchild), _dptr(F), _dptr(T)),
               "pr_mlp_features")
        return F, T

    def mlp_warm_start(self, nodes, params, Bparent):
        """(B0, choice, gaps): starting points for child nodes, the FP64 gap
        deciding between the parent solution (choice 0), prox(beta_parent)
        (1) and, with params, the network's candidate (2); gaps (m, 3) in that
        order."""
        import torch
        m = len(nodes)
        dev = self.X.device
        arr = (PrNode * m)(*[nd.c() for nd in nodes])
        Bparent = Bparent.to(device=dev, dtype=torch.float64).contiguous()
        B0 = torch.empty_like(Bparent)
        choice = (ctypes.c_int32 * max(m, 1))()
        gaps = (ctypes.c_double * max(3 * m, 1))()
        _check(load().pr_mlp_warm_start(self.h, arr, m, _dptr(None if params is None else params.contiguous()),
                                        _dptr(Bparent), _dptr(B0), choice, gaps), "pr_mlp_warm_start")
        return B0, np.array(choice[:m], dtype=np.int32), np.array(gaps[:3 * m]).reshape(m, 3)

    def dual_bound(self, node, zeta=None, beta=None):
        lb = ctypes.c_double()
        ph = ctypes.c_double(float("nan"))
        nd = node.c()
        _check(load().pr_dual_bound(self.h, ctypes.byref(nd), _dptr(zeta), _dptr(beta), ctypes.byref(lb),
                                    ctypes.byref(ph)), "pr_dual_bound")
        return lb.value, ph.value

    def gemv(self, b):
        import torch
        u = torch.empty(self.n, dtype=torch.float64, device=self.X.device)
        _check(load().pr_gemv(self.h, _dptr(b.contiguous()), _dptr(u)), "pr_gemv")
        return u

    def gemv_t(self, r):
        import torch
        h = torch.empty(self.p, dtype=torch.float64, device=self.X.device)
        _check(load().pr_gemv_t(self.h, _dptr(r.contiguous()), _dptr(h)), "pr_gemv_t")
        return h

    def gemv_t2(self, r1, r2):
        import torch
        h1 = torch.empty(self.p, dtype=torch.float64, device=self.X.device)
        h2 = torch.empty(self.p, dtype=torch.float64, device=self.X.device)
        _check(load().pr_gemv_t2(self.h, _dptr(r1.contiguous()), _dptr(r2.contiguous()), _dptr(h1), _dptr(h2)),
               "pr_gemv_t2")
        return h1, h2

    def time_gemv(self, b, reps=20):
        import torch
        u = torch.empty(self.n, dtype=torch.float64, device=self.X.device)
        ms = ctypes.c_double()
        _check(load().pr_time_gemv(self.h, _dptr(b.contiguous()), _dptr(u), int(reps), ctypes.byref(ms)),
               "pr_time_gemv")
        return ms.value

    def time_gemv_t(self, r, reps=20):
        import torch
        h = torch.empty(self.p, dtype=torch.float64, device=self.X.device)
        ms = ctypes.c_double()
        _check(load().pr_time_gemv_t(self.h, _dptr(r.contiguous()), _dptr(h), int(reps), ctypes.byref(ms)),
               "pr_time_gemv_t")
        return ms.value


def prox(v, rho, k, M, status):
    """prox_{rho g_N}(v) on the device (v: CUDA float64, status: CUDA int8)."""
    import torch
    out = torch.empty_like(v)
    _check(load().pr_prox(_stream_ptr(), _dptr(v.contiguous()), v.numel(), float(rho), int(k), float(M),
                          _dptr(status.contiguous()), _dptr(out)), "pr_prox")
    return out


def prox_noalloc(v, rho, k, M, status, out=None):
    """prox_{rho g_N}(v) through pr_prox_noalloc (no allocation inside the
    library; `out`, a CUDA float64 tensor like v, is allocated here if not
    given)."""
    import torch
    if out is None:
        out = torch.empty_like(v)
    _check(load().pr_prox_noalloc(_stream_ptr(), _dptr(v.contiguous()), v.numel(), float(rho), int(k), float(M),
                                  _dptr(status.contiguous()), _dptr(out)), "pr_prox_noalloc")
    return out


def time_prox(v, rho, k, M, status, reps=20):
    """(prox output, ms per prox launch, ms per g_N launch) on the device."""
    import torch
    out = torch.empty_like(v)
    a = ctypes.c_double()
    b = ctypes.c_double()
    _check(load().pr_time_prox(_stream_ptr(), _dptr(v.contiguous()), v.numel(), float(rho), int(k), float(M),
                               _dptr(status.contiguous()), _dptr(out), int(reps), ctypes.byref(a), ctypes.byref(b)),
           "pr_time_prox")
    return out, a.value, b.value


def time_read(buf, blocks, unroll=1, reps=20):
    """ms per plain streaming read of the CUDA tensor `buf` (pr_time_read,
    on the current stream)."""
    ms = ctypes.c_double()
    _check(load().pr_time_read(_dptr(buf), buf.numel() * buf.element_size(), int(blocks), int(unroll), int(reps),
                               _stream_ptr(), ctypes.byref(ms)), "pr_time_read")
    return ms.value


def gemm(A, B, KS=1):
    """C[z] = B[:, split z] @ A[:, split z]^T for a bfloat16 CUDA tensor A
    (Mc x K) and a float64 CUDA tensor B (Nr x K), FP64 MFMA; returns
    (KS, Nr, Mc) float64."""
    import torch
    if A.dtype != torch.bfloat16 or B.dtype != torch.float64 or A.stride(1) != 1 or B.stride(1) != 1:
        raise ValueError("gemm: A bfloat16 and B float64, both row-major")
    Mc, K = A.shape
    Nr = B.shape[0]
    C = torch.empty((KS, Nr, Mc), dtype=torch.float64, device=A.device)
    _check(load().pr_gemm(_stream_ptr(), _dptr(A), A.stride(0), _dptr(B), B.stride(0), _dptr(C), Mc, Nr, K, int(KS)),
           "pr_gemm")
    return C


def mlp_forward(params, F):
    """Network output (rows,) float32 for feature rows F (rows, 8) bfloat16."""
    import torch
    out = torch.empty(F.shape[0], dtype=torch.float32, device=F.device)
    _check(load().pr_mlp_forward(_stream_ptr(), _dptr(params), _dptr(F.contiguous()), F.shape[0], _dptr(out)),
           "pr_mlp_forward")
    return out


def mlp_workspace(rows):
    return int(load().pr_mlp_workspace(int(rows)))


def mlp_grad(params, F, T, work=None, grad=None):
    """(gradient (4801,), loss) of the mean squared error; work / grad may be
    preallocated float32 device tensors of mlp_workspace(rows) / 4802 entries."""
    import torch
    rows = F.shape[0]
    if work is None:
        work = torch.empty(mlp_workspace(rows), dtype=torch.float32, device=F.device)
    if grad is None:
        grad = torch.empty(MLP_NPARAM + 1, dtype=torch.float32, device=F.device)
    _check(load().pr_mlp_grad(_stream_ptr(), _dptr(params), _dptr(F), _dptr(T), rows, _dptr(work), _dptr(grad)),
           "pr_mlp_grad")
    return grad


def mlp_adam(params, grad, m1, m2, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on params (float32 device) from grad[:4801]."""
    _check(load().pr_mlp_adam(_stream_ptr(), _dptr(params), _dptr(grad), _dptr(m1), _dptr(m2), int(step),
                              float(lr), float(beta1), float(beta2), float(eps)), "pr_mlp_adam")


def regularizer(beta, alpha, k, M, status):
    """(g_N(beta), g_N*(alpha)) computed on the device; either input may be None."""
    g = ctypes.c_double(float("nan"))
    gs = ctypes.c_double(float("nan"))
    p = (beta if beta is not None else alpha).numel()
    _check(load().pr_regularizer(_stream_ptr(), _dptr(beta), _dptr(alpha), p, int(k), float(M),
                                 _dptr(status.contiguous()),
                                 ctypes.byref(g) if beta is not None else None,
                                 ctypes.byref(gs) if alpha is not None else None), "pr_regularizer")
    return (g.value if beta is not None else None, gs.value if alpha is not None else None)


E3 = math.exp(3.0)
