"""Learned warm start for child nodes: training data from a seeded random
branching process, training of the per-coordinate network, and its
evaluation against the parent warm start.

Control flow only: every arithmetic step (node solves, feature rows, network
forward and backward, Adam, the FP64 gap that accepts or rejects a proposal)
runs in libpr's kernels; torch holds device memory and gathers rows.

Branching process: a pool of solved nodes starts at the root; each round draws
m parents uniformly from the pool, branches each on a uniformly random free
coordinate, fixed to one or to zero by a fair coin (to zero when the parent
already fixes k coordinates to one), and solves the m children together with
the parents' solutions as starting points.  Each child gives one training pair
(parent solution, child solution), i.e. p feature rows with targets
beta_child - beta_parent, and joins the pool.
"""
import time

import numpy as np

from ._binding import Node, FREE, CONVERGED, MLP_NFEAT, MLP_NPARAM, mlp_grad, mlp_adam, mlp_workspace

H = 64


def init_params(seed, device):
    """He-uniform weights (bound sqrt(6 / fan_in)), output layer scaled by 0.1,
    zero biases; float32 on `device`."""
    import torch
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, MLP_NFEAT)) * np.sqrt(6.0 / MLP_NFEAT)
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    w3 = rng.uniform(-1, 1, H) * np.sqrt(6.0 / H) * 0.1
    P = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, [0.0]])
    assert P.size == MLP_NPARAM
    return torch.tensor(P, dtype=torch.float32, device=device)


def random_children(parents, p, rng):
    """One child per parent, branched on a uniformly random free coordinate."""
    out = []
    for nd in parents:
        free = np.flatnonzero(nd.status(p) == FREE)
        j = int(free[rng.integers(free.size)])
        if rng.random() < 0.5 and nd.J1.size < nd.k:
            out.append(Node(nd.k, nd.lambda2, nd.M, J0=nd.J0, J1=np.append(nd.J1, j)))
        else:
            out.append(Node(nd.k, nd.lambda2, nd.M, J0=np.append(nd.J0, j), J1=nd.J1))
    return out


class BranchingPool:
    """Solved nodes of the branching process; their solutions stay on the device."""

    def __init__(self, ctx, root, capacity, **opts):
        import torch
        self.ctx = ctx
        self.p = ctx.p
        self.opts = opts
        self.B = torch.empty((capacity, self.p), dtype=torch.float64, device=ctx.X.device)
        res, B = ctx.solve_batch([root], **opts)
        if res[0]["status"] != CONVERGED:
            raise RuntimeError(f"root solve did not converge: {res[0]}")
        self.B[0].copy_(B[0])
        self.nodes = [root]

    def grow(self, m, rng, keep=True):
        """Branch m uniformly drawn parents once each and solve the children;
        returns (children, parent solutions (m, p), child solutions (m, p), results)."""
        import torch
        idx = rng.integers(0, len(self.nodes), m)
        children = random_children([self.nodes[i] for i in idx], self.p, rng)
        Bp = self.B[torch.as_tensor(idx, device=self.B.device)]
        res, Bc = self.ctx.solve_batch(children, B0=Bp, **self.opts)
        if keep:
            n0 = len(self.nodes)
            take = min(m, self.B.shape[0] - n0)
            if take > 0:
                self.B[n0:n0 + take].copy_(Bc[:take])
                self.nodes.extend(children[:take])
        return children, Bp, Bc, res


def generate_pairs(pool, n_pairs, batch, rng, progress=None):
    """Feature rows F (n_pairs * p, 8) bfloat16 and targets T (n_pairs * p,)
    float32 from n_pairs children of the branching process."""
    import torch
    p = pool.p
    dev = pool.B.device
    F = torch.empty((n_pairs * p, MLP_NFEAT), dtype=torch.bfloat16, device=dev)
    T = torch.empty(n_pairs * p, dtype=torch.float32, device=dev)
    done = 0
    iters = []
    while done < n_pairs:
        m = min(batch, n_pairs - done)
        children, Bp, Bc, res = pool.grow(m, rng)
        f, t = pool.ctx.mlp_features(children, Bp, Bc)
        F[done * p:(done + m) * p].copy_(f)
        T[done * p:(done + m) * p].copy_(t)
        iters.extend(r["iters"] for r in res)
        done += m
        if progress:
            progress(done, n_pairs)
    return F, T, np.array(iters)


def train(params, F, T, epochs, batch_rows, lr, seed, progress=None):
    """Adam on the mean squared error over minibatches of batch_rows
    consecutive rows, in a fresh random order every epoch.  Returns the mean
    minibatch loss of every epoch."""
    import torch
    rows = F.shape[0]
    nb = max(1, rows // batch_rows)
    dev = F.device
    work = torch.empty(mlp_workspace(batch_rows), dtype=torch.float32, device=dev)
    grad = torch.empty(MLP_NPARAM + 1, dtype=torch.float32, device=dev)
    m1 = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev)
    m2 = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev)
    hist = torch.empty(nb, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    losses = []
    step = 0
    for ep in range(epochs):
        for q, b in enumerate(rng.permutation(nb)):
            r0 = int(b) * batch_rows
            r1 = rows if b == nb - 1 else r0 + batch_rows
            if r1 - r0 != batch_rows:
                w = torch.empty(mlp_workspace(r1 - r0), dtype=torch.float32, device=dev)
            else:
                w = work
            mlp_grad(params, F[r0:r1], T[r0:r1], w, grad)
            step += 1
            mlp_adam(params, grad, m1, m2, step, lr=lr)
            hist[q].copy_(grad[MLP_NPARAM])
        losses.append(float(np.mean(hist.cpu().numpy().astype(np.float64))))
        if progress:
            progress(ep, losses[-1])
    return losses


def _solve_chunks(ctx, children, B0, **opts):
    res = []
    for a in range(0, len(children), ctx.max_batch):
        r, _ = ctx.solve_batch(children[a:a + ctx.max_batch], B0=B0[a:a + ctx.max_batch], want_beta=False, **opts)
        res.extend(r)
    return res


def evaluate(ctx, params, children, Bp, **opts):
    """Iterations and wall time to the FP64 gap tolerance from three starts:
    the parent solutions, the judged start without the network (the smaller
    FP64 gap of the parent and prox(beta_parent); pr_mlp_warm_start with no
    parameters) and the judged start with it (the smallest gap of those two
    and prox(beta_parent + output)).  Times of the judged starts include
    building them."""
    import torch

    def run(make_start):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B0, choice, gaps = make_start()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = _solve_chunks(ctx, children, B0, **opts)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return res, t1 - t0, t2 - t1, choice, gaps

    rp, _, sp, _, _ = run(lambda: (Bp, None, None))
    ra, wa, sa, ca, ga = run(lambda: ctx.mlp_warm_start(children, None, Bp))
    rm, wm, sm, cm, gm = run(lambda: ctx.mlp_warm_start(children, params, Bp))
    ip = np.array([r["iters"] for r in rp])
    ia = np.array([r["iters"] for r in ra])
    im = np.array([r["iters"] for r in rm])
    ok = all(r["status"] == CONVERGED for rr in (rp, ra, rm) for r in rr)

    def bound_diff(x):
        return float(max(abs(a["lower_bound"] - b["lower_bound"]) / abs(a["primal"]) for a, b in zip(rp, x)))

    return {"nodes": len(children), "all_converged": ok,
            "parent_iters_mean": float(ip.mean()), "parent_iters_median": float(np.median(ip)),
            "prox_parent_iters_mean": float(ia.mean()), "prox_parent_iters_median": float(np.median(ia)),
            "learned_iters_mean": float(im.mean()), "learned_iters_median": float(np.median(im)),
            "parent_solve_s": sp,
            "prox_parent_start_s": wa, "prox_parent_solve_s": sa, "prox_parent_total_s": wa + sa,
            "learned_start_s": wm, "learned_solve_s": sm, "learned_total_s": wm + sm,
            "prox_parent_start_kept": float(np.mean(ca == 1)), "network_start_kept": float(np.mean(cm == 2)),
            "parent_gap_median": float(np.median(gm[:, 0])),
            "prox_parent_start_gap_median": float(np.median(np.min(ga[:, :2], axis=1))),
            "learned_start_gap_median": float(np.median(np.min(gm, axis=1))),
            "max_rel_bound_difference": max(bound_diff(ra), bound_diff(rm)),
            "iters_parent": ip, "iters_prox_parent": ia, "iters_learned": im, "choice": cm, "gaps": gm}
