"""Learned warm start on the GPU: the network's forward pass, gradient and
Adam step against the FP64 oracle, the feature rows against the oracle's
features, the FP64-gap judge of pr_mlp_warm_start, and what a trained network
gains over the parent warm start on a small branching process.

Tolerances.  The kernels round the weights, the features' products and the
hidden activations to BF16 (relative error <= 2^-8 each) and accumulate in
FP32; the oracle computes in FP64 from the FP32 master weights.  The forward
bound below propagates those roundings through absolute values of the
oracle's own layers; gradients are products of at most four rounded factors,
so each entry is within about 4 * 2^-8 relative of its terms, checked as a
2.5% bound on each parameter block's norm."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from workloads import make_instance

pytestmark = pytest.mark.gpu

U = 2.0 ** -8      # BF16 unit roundoff (8-bit significand)


def _pr():
    import paper_2603_01306_amd as pr
    return pr


def _bf16(a):
    """Round float64 values to the nearest BF16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((f + 0x7FFF + ((f >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _rand_params(seed, bf16_weights=True):
    """FP32 master values; with bf16_weights the matrix weights W1, W2 are
    BF16 numbers, so the kernels' weight rounding is exact and a ReLU mask can
    only differ where a pre-activation is within FP32 rounding of zero."""
    rng = np.random.default_rng(seed)
    P = omlp.init_params(seed)
    P[omlp.OFF_B1:omlp.OFF_W2] = rng.normal(0, 0.3, omlp.H)
    P[omlp.OFF_B2:omlp.OFF_W3] = rng.normal(0, 0.3, omlp.H)
    P[omlp.OFF_W3:omlp.OFF_B3] *= 10.0
    P[omlp.OFF_B3] = 0.1
    if bf16_weights:
        P[omlp.OFF_W1:omlp.OFF_B1] = _bf16(P[omlp.OFF_W1:omlp.OFF_B1])
        P[omlp.OFF_W2:omlp.OFF_B2] = _bf16(P[omlp.OFF_W2:omlp.OFF_B2])
    return P.astype(np.float32).astype(np.float64)


def _rand_rows(seed, rows):
    rng = np.random.default_rng(seed)
    F = _bf16(rng.normal(0, 1, (rows, omlp.NF)))
    T = rng.normal(0, 1, rows).astype(np.float32).astype(np.float64)
    return F, T


def _dev(a, dt):
    import torch
    return torch.tensor(a, dtype=dt, device="cuda")


def _forward_bound(P, F):
    """First-order bound on |out_gpu - out_oracle| from BF16 rounding of W1,
    W2, a1 and the FP32 sums, propagated through absolute values (x2 margin)."""
    W1, b1, W2, b2, w3, b3 = omlp.unpack(P)
    A = np.abs(F) @ np.abs(W1).T
    z1 = F @ W1.T + b1
    e1 = U * A + 1e-6 * (A + np.abs(b1))
    a1 = np.maximum(z1, 0)
    e1 = e1 + U * np.abs(a1)
    e2 = e1 @ np.abs(W2).T + U * (np.abs(a1) @ np.abs(W2).T) + 1e-6 * (np.abs(a1) @ np.abs(W2).T + np.abs(b2))
    return 2.0 * (e2 @ np.abs(w3)) + 1e-6


@pytest.mark.parametrize("rows", [1, 31, 3000, 131109])
def test_forward_matches_oracle(dev, rows):
    import torch
    pr = _pr()
    P = _rand_params(rows, bf16_weights=rows % 2 == 1)
    F, _ = _rand_rows(rows + 1, rows)
    out = pr.mlp_forward(_dev(P, torch.float32), _dev(F, torch.float32).to(torch.bfloat16)).cpu().numpy()
    ref = omlp.forward(P, F)
    assert np.all(np.abs(out - ref) <= _forward_bound(P, F))


@pytest.mark.parametrize("rows", [37, 5000, 131109])
def test_gradient_matches_oracle(dev, rows):
    """131109 rows take several row chunks per workgroup and a ragged tail."""
    import torch
    pr = _pr()
    P = _rand_params(7 + rows)
    F, T = _rand_rows(9 + rows, rows)
    g = pr.mlp_grad(_dev(P, torch.float32), _dev(F, torch.float32).to(torch.bfloat16),
                    _dev(T, torch.float32)).cpu().numpy().astype(np.float64)
    loss, ref = omlp.loss_grad(P, F, T)
    assert abs(g[-1] - loss) <= 0.02 * loss
    blocks = [(omlp.OFF_W1, omlp.OFF_B1), (omlp.OFF_B1, omlp.OFF_W2), (omlp.OFF_W2, omlp.OFF_B2),
              (omlp.OFF_B2, omlp.OFF_W3), (omlp.OFF_W3, omlp.OFF_B3), (omlp.OFF_B3, omlp.NPARAM)]
    for a, b in blocks:
        err = np.linalg.norm(g[a:b] - ref[a:b])
        assert err <= 0.025 * np.linalg.norm(ref[a:b]) + 1e-7, (a, b, err, np.linalg.norm(ref[a:b]))


def _grad_error_bound(P, F, T):
    """Per-parameter bound on |g_gpu - g_oracle(P_bf16)| where P_bf16 rounds
    W1, W2 to BF16 as the kernels do.  Errors are propagated through absolute
    values of the oracle's own layers: FP32 accumulation (1e-6 of the absolute
    sum), BF16 rounding (U) of a1 and of dz2, dz1 where they enter an MFMA
    product, and every ReLU mask whose pre-activation is within its own error
    bound of zero counted as fully uncertain.  A factor 2 covers second-order
    terms."""
    W1, b1, W2, b2, w3, b3 = omlp.unpack(P)
    N = F.shape[0]
    aF, aW1, aW2, aw3 = np.abs(F), np.abs(W1), np.abs(W2), np.abs(w3)
    eps32 = 1e-6
    z1 = F @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    Ez1 = eps32 * (aF @ aW1.T + np.abs(b1))
    Ea1 = Ez1 + U * a1
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    Ez2 = Ea1 @ aW2.T + eps32 * (a1 @ aW2.T + np.abs(b2))
    Ea2 = Ez2 + U * a2
    out = a2 @ w3 + b3
    Eout = Ea2 @ aw3 + eps32 * (a2 @ aw3 + abs(b3))
    dout = 2.0 * (out - T) / N
    Edout = 2.0 * Eout / N
    u1, u2 = np.abs(z1) <= Ez1, np.abs(z2) <= Ez2          # masks that may flip
    dz2 = np.outer(dout, w3) * (z2 > 0)
    Edz2 = np.outer(Edout, aw3) + U * np.abs(dz2) + u2 * np.abs(np.outer(dout, w3))
    dz1 = (dz2 @ W2) * (z1 > 0)
    Edz1 = (Edz2 @ aW2 + U * (np.abs(dz2) @ aW2)) * ((z1 > 0) | u1) + u1 * (np.abs(dz2) @ aW2)
    gW3 = Edout @ a2 + np.abs(dout) @ Ea2 + eps32 * (np.abs(dout) @ a2)
    gB3 = np.sum(Edout) + eps32 * np.sum(np.abs(dout))
    gW2 = Edz2.T @ a1 + np.abs(dz2).T @ Ea1 + eps32 * (np.abs(dz2).T @ a1)
    gB2 = Edz2.sum(axis=0) + eps32 * np.abs(dz2).sum(axis=0)
    gW1 = Edz1.T @ aF + eps32 * (np.abs(dz1).T @ aF)
    gB1 = Edz1.sum(axis=0) + eps32 * np.abs(dz1).sum(axis=0)
    return 2.0 * omlp.pack(gW1, gB1, gW2, gB2, gW3, gB3) + 1e-9


@pytest.mark.parametrize("rows", [37, 5000, 131109])
def test_gradient_with_fp32_master_weights(dev, rows):
    """General FP32 master weights (training's case, not BF16-exact): each
    gradient entry against the oracle evaluated at the BF16-rounded weights
    the kernels use, within a bound derived per entry from the arithmetic."""
    import torch
    pr = _pr()
    P = _rand_params(11 + rows, bf16_weights=False)
    F, T = _rand_rows(13 + rows, rows)
    Pb = P.copy()
    Pb[omlp.OFF_W1:omlp.OFF_B1] = _bf16(P[omlp.OFF_W1:omlp.OFF_B1])
    Pb[omlp.OFF_W2:omlp.OFF_B2] = _bf16(P[omlp.OFF_W2:omlp.OFF_B2])
    assert np.any(Pb != P)
    g = pr.mlp_grad(_dev(P, torch.float32), _dev(F, torch.float32).to(torch.bfloat16),
                    _dev(T, torch.float32)).cpu().numpy().astype(np.float64)
    loss, ref = omlp.loss_grad(Pb, F, T)
    bound = _grad_error_bound(Pb, F, T)
    err = np.abs(g[:-1] - ref)
    worst = int(np.argmax(err / bound))
    print(f"rows={rows} max err/bound={err[worst] / bound[worst]:.3f} at {worst}, "
          f"median bound/|g|={np.median(bound / (np.abs(ref) + 1e-30)):.3g}", flush=True)
    assert np.all(err <= bound), (worst, err[worst], bound[worst], ref[worst])
    assert abs(g[-1] - loss) <= 0.02 * loss
    # the entry bounds grow where a gradient sums terms of both signs; each
    # parameter block as a whole stays within a few BF16 roundings
    blocks = [(omlp.OFF_W1, omlp.OFF_B1), (omlp.OFF_B1, omlp.OFF_W2), (omlp.OFF_W2, omlp.OFF_B2),
              (omlp.OFF_B2, omlp.OFF_W3), (omlp.OFF_W3, omlp.OFF_B3), (omlp.OFF_B3, omlp.NPARAM)]
    for a, b in blocks:
        rel = np.linalg.norm(g[a:b] - ref[a:b]) / (np.linalg.norm(ref[a:b]) + 1e-30)
        print(f"  block {a}:{b} relative error {rel:.2e}", flush=True)
        assert rel <= 0.025


def test_gradient_is_deterministic(dev):
    import torch
    pr = _pr()
    P = _dev(_rand_params(3), torch.float32)
    F, T = _rand_rows(4, 70000)
    Fd, Td = _dev(F, torch.float32).to(torch.bfloat16), _dev(T, torch.float32)
    assert torch.equal(pr.mlp_grad(P, Fd, Td), pr.mlp_grad(P, Fd, Td))


def test_adam_matches_oracle(dev):
    import torch
    pr = _pr()
    rng = np.random.default_rng(5)
    P = rng.normal(size=omlp.NPARAM).astype(np.float32).astype(np.float64)
    Pd = _dev(P, torch.float32)
    m1 = torch.zeros(omlp.NPARAM, dtype=torch.float32, device="cuda")
    m2 = torch.zeros_like(m1)
    m, v = np.zeros(omlp.NPARAM), np.zeros(omlp.NPARAM)
    for step in range(1, 6):
        g = rng.normal(size=omlp.NPARAM + 1).astype(np.float32).astype(np.float64)
        pr.mlp_adam(Pd, _dev(g, torch.float32), m1, m2, step, lr=0.01)
        P, m, v = omlp.adam(P, g[:-1], m, v, step, lr=0.01)
    assert np.allclose(Pd.cpu().numpy(), P, rtol=1e-6, atol=1e-6)


@pytest.fixture(scope="module")
def inst_ctx(dev):
    import torch
    pr = _pr()
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=0, seed=31, storage="bf16")
    X = torch.from_numpy(inst.Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
    ctx = pr.Context(X, torch.from_numpy(inst.y).to(dev), 0, max_batch=64)
    yield inst, ctx
    ctx.close()


def test_features_match_oracle(inst_ctx):
    import torch
    pr = _pr()
    inst, ctx = inst_ctx
    rng = np.random.default_rng(11)
    nodes = [pr.Node(8, 0.2, 2.0, J0=[3, 40], J1=[7]), pr.Node(8, 0.2, 2.0), pr.Node(5, 0.5, 2.0, J1=[1, 2])]
    Bp = np.zeros((3, inst.p))
    for i in range(3):
        nz = rng.choice(inst.p, 12, replace=False)
        Bp[i, nz] = rng.normal(size=12)
    Bp[1, 5] = Bp[1, 9] = 0.75                    # tied magnitudes
    Bc = Bp + rng.normal(0, 0.01, Bp.shape)
    F, T = ctx.mlp_features(nodes, torch.tensor(Bp, device="cuda"), torch.tensor(Bc, device="cuda"))
    F = F.float().cpu().numpy().astype(np.float64).reshape(3, inst.p, 8)
    T = T.cpu().numpy().reshape(3, inst.p)
    X = inst.X64().T                  # (n, p)
    for i, nd in enumerate(nodes):
        st = nd.status(inst.p)
        w = oracle.rmatvec(inst.Xcm, 2.0 * (inst.y - X @ Bp[i]))      # X^T zeta at the parent
        ref = omlp.features(Bp[i], w, st, nd.lambda2, nd.k)
        # one BF16 rounding of FP64 values (the GPU rounds through FP32)
        assert np.all(np.abs(F[i] - _bf16(ref)) <= 2 * U * np.abs(ref) + 1e-30)
        assert np.array_equal(T[i], (Bc[i] - Bp[i]).astype(np.float32))


@pytest.mark.parametrize("batched", [True, False])
@pytest.mark.parametrize("with_net", [True, False])
def test_warm_start_judge(inst_ctx, dev, batched, with_net):
    """Every reported gap is the oracle's FP64 gap of its candidate (the parent,
    prox(beta_parent) -- exactly the oracle's prox_{rho g_N} with rho =
    2 lambda2 / L -- and, with a network, its proposal), and the start kept is
    the candidate with the smallest gap; the batched evaluation (all children
    at once) and the one-at-a-time path alike."""
    import torch
    pr = _pr()
    inst, bctx = inst_ctx
    from paper_2603_01306_amd import learned
    if batched:
        ctx = bctx
    else:
        X = torch.from_numpy(inst.Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
        ctx = pr.Context(X, torch.from_numpy(inst.y).to(dev), 0, max_batch=1)
    rng = np.random.default_rng(2)
    root = pr.Node(8, 0.2, 2.0)
    res, Br = ctx.solve_batch([root], rel_gap_tol=1e-8)
    children = learned.random_children([root] * 6, inst.p, rng)
    children.append(pr.Node(2, 0.2, 2.0, J1=[1, 2, 3]))       # infeasible: keeps the parent
    Bp = Br.repeat(len(children), 1)
    params = learned.init_params(0, "cuda") if with_net else None
    B0, choice, gaps = ctx.mlp_warm_start(children, params, Bp)
    B0 = B0.cpu().numpy()
    L = 1.01 * 2.0 * ctx.norm2()
    X = inst.X64().T

    def gap(st, b):
        ph = oracle.primal(inst.Xcm, inst.y, b, 0, 0.2, 2.0, 8, status=st)
        if not math.isfinite(ph):
            return math.inf, ph
        zeta = 2.0 * (inst.y - X @ b)
        return ph - oracle.dual(inst.Xcm, inst.y, zeta, 0, 0.2, 2.0, 8, status=st), ph

    for i, nd in enumerate(children):
        st = nd.status(inst.p)
        par = Bp[i].cpu().numpy()
        if i == len(children) - 1:
            assert choice[i] == 0 and np.array_equal(B0[i], par) and np.all(np.isinf(gaps[i]))
            continue
        assert choice[i] == int(np.argmin(gaps[i]))
        if not with_net:
            assert math.isinf(gaps[i, 2])
        gp, php = gap(st, par)
        assert (math.isinf(gp) and math.isinf(gaps[i, 0])) or abs(gp - gaps[i, 0]) <= 1e-9 * abs(php)
        pp = oracle.prox_g(par, 2.0 * 0.2 / L, 8, 2.0, st)
        ga, pha = gap(st, pp)
        assert abs(ga - gaps[i, 1]) <= 1e-9 * abs(pha)
        if choice[i] == 0:
            assert np.array_equal(B0[i], par)
        elif choice[i] == 1:
            assert np.max(np.abs(B0[i] - pp)) <= 1e-12 * max(1.0, np.max(np.abs(pp)))
        else:
            gn, phn = gap(st, B0[i])
            assert abs(gn - gaps[i, 2]) <= 1e-9 * abs(phn)
    assert np.sum(choice[:-1] > 0) >= 1
    if not batched:
        ctx.close()


def test_training_gains_over_parent_start(inst_ctx):
    """Train on children of a small branching process; on held-out children
    the network predicts the child solutions better than the parent solution
    does (lower mean squared error of the warm start), and solving from the
    judged starts reaches the same bounds."""
    import torch
    pr = _pr()
    from paper_2603_01306_amd import learned
    inst, ctx = inst_ctx
    rng = np.random.default_rng(4)
    pool = learned.BranchingPool(ctx, pr.Node(8, 0.2, 2.0), capacity=1200, rel_gap_tol=1e-7)
    F, T, it = learned.generate_pairs(pool, 640, 64, rng)
    params = learned.init_params(1, "cuda")
    losses = learned.train(params, F, T, epochs=12, batch_rows=8192, lr=2e-3, seed=3)
    print("losses", [round(x, 6) for x in losses], flush=True)
    assert losses[-1] < losses[0]
    children, Bp, Bc, _ = pool.grow(64, rng, keep=False)
    Fh, Th = ctx.mlp_features(children, Bp, Bc)
    out = pr.mlp_forward(params, Fh)
    mse_net = float(np.mean((out.cpu().numpy().astype(np.float64) - Th.cpu().numpy()) ** 2))
    mse_par = float(np.mean(Th.cpu().numpy().astype(np.float64) ** 2))
    print("held-out mse: network", mse_net, "parent", mse_par, flush=True)
    assert mse_net < mse_par
    ev = learned.evaluate(ctx, params, children, Bp, rel_gap_tol=1e-7)
    print({k: v for k, v in ev.items() if not isinstance(v, np.ndarray)}, flush=True)
    assert ev["all_converged"] and ev["max_rel_bound_difference"] <= 2e-7
    # what the network adds over the same judged start without it: its
    # candidate joins the judged ones, so the start gap can only fall; the
    # held-out iterations of the three starts are reported (the gain is small,
    # and on this branching process the network's candidate is rarely kept)
    print("iterations: parent", ev["parent_iters_mean"], "prox(parent)", ev["prox_parent_iters_mean"],
          "network", ev["learned_iters_mean"], "network kept", ev["network_start_kept"], flush=True)
    assert ev["learned_start_gap_median"] <= ev["prox_parent_start_gap_median"]
    assert ev["prox_parent_start_gap_median"] <= ev["parent_gap_median"]
