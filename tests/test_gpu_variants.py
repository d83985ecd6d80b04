"""AC-FGM (with and without the duality-gap restart) and the LASSO solves with
the gap restart on the GPU, through the C ABI, against the oracle: the
per-evaluation (Phi, Psi) traces, iteration / restart / line-search counts,
and at full size the certificates recomputed by the oracle."""
import math

import numpy as np
import pytest

import oracle
from workloads import make_instance, config_instance

pytestmark = pytest.mark.gpu


def _ctx(dev, inst):
    import torch
    import paper_2603_01306_amd as pr
    return pr.Context(torch.from_numpy(inst.Xcm).to(dev), torch.from_numpy(inst.y).to(dev), inst.loss)


def _trace(dev, its):
    import torch
    return torch.full((2 * (its + 1),), float("nan"), dtype=torch.float64, device=dev)


@pytest.mark.parametrize("loss,storage,restart", [(0, "f64", True), (0, "f32", False), (1, "f64", True),
                                                  (1, "f32", False)])
def test_acfgm_trace_matches_oracle(dev, loss, storage, restart):
    import paper_2603_01306_amd as pr
    inst = make_instance(n=512, p=200, corr=0.6, k_true=6, snr=5.0, loss=loss, seed=50 + loss, storage=storage)
    ctx = _ctx(dev, inst)
    node = pr.Node(6, 0.4, 2.0, J0=[3, 17], J1=[8])
    st = node.status(inst.p)
    L = (2.0 if loss == 0 else 0.25) * float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max()) * 1.01
    L0, its = L / 40.0, 300
    tr = _trace(dev, its)
    method = pr.ACFGM_GAP if restart else pr.ACFGM
    r = ctx.solve(node, want_zeta=True, rel_gap_tol=1e-9, max_iter=its, L0=L0, acfgm_b=0.1, acfgm_c=2.0,
                  method=method, eta=math.e, trace=tr)
    ref = oracle.solve_acfgm(inst.Xcm, inst.y, loss, 0.4, 2.0, 6, status=st, L0=L0, c=2.0, b=0.1, restart=restart,
                             tol=1e-9, eta=math.e, max_iter=its, trace_cap=its + 1)
    print({k: v for k, v in r.items() if k not in ("beta", "zeta")}, ref["iters"], ref["restarts"], ref["rejected"],
          flush=True)
    assert r["iters"] == ref["iters"] and r["restarts"] == ref["restarts"] and r["trials"] == ref["rejected"]
    assert r["trials"] >= 1 and r["L"] == pytest.approx(ref["L1"], rel=1e-15)
    t = tr.cpu().numpy().reshape(-1, 2)[: r["iters"] + 1]
    scale = abs(ref["ub"])
    np.testing.assert_allclose(t[:, 0], ref["phi_trace"], rtol=0, atol=1e-10 * scale)
    np.testing.assert_allclose(t[:, 1], ref["phi_trace"] - ref["trace"], rtol=0, atol=1e-10 * scale)
    assert abs(r["lower_bound"] - ref["lb"]) <= 1e-10 * scale and abs(r["primal"] - ref["ub"]) <= 1e-10 * scale
    psi = oracle.dual(inst.Xcm, inst.y, r["zeta"].cpu().numpy(), loss, 0.4, 2.0, 6, status=st)
    assert abs(psi - r["lower_bound"]) <= 1e-12 * scale
    phi = oracle.primal(inst.Xcm, inst.y, r["beta"].cpu().numpy(), loss, 0.4, 2.0, 6, status=st)
    assert abs(phi - r["primal"]) <= 1e-12 * scale
    ctx.close()


def test_acfgm_gap_restart_converges_on_the_full_size_root(dev):
    """n = 16384, p = 8192 FP32 least-squares root with AC-FGM + gap restart to
    1e-6: the certificate (zeta, beta) recomputed over the stored X."""
    import paper_2603_01306_amd as pr
    inst = config_instance("ls_root_n16384_p8192_f32")
    ctx = _ctx(dev, inst)
    r = ctx.solve(pr.Node(20, 0.1, 2.0), want_zeta=True, method=pr.ACFGM_GAP, max_iter=20000)
    print({k: v for k, v in r.items() if k not in ("beta", "zeta")}, flush=True)
    assert r["status"] == pr.CONVERGED and r["restarts"] >= 3
    psi = oracle.dual(inst.Xcm, inst.y, r["zeta"].cpu().numpy(), 0, 0.1, 2.0, 20)
    phi = oracle.primal(inst.Xcm, inst.y, r["beta"].cpu().numpy(), 0, 0.1, 2.0, 20)
    assert abs(psi - r["lower_bound"]) <= 1e-10 * abs(psi)
    assert abs(phi - r["primal"]) <= 1e-10 * abs(phi)
    assert 0.0 <= (phi - psi) / abs(phi) <= 1e-6
    ctx.close()


def _lam(inst, kind, frac):
    X = inst.X64().T
    if kind == oracle.L1_REG:
        return frac * 2.0 * float(np.max(np.abs(X.T @ inst.y)))   # a fraction of the smallest lam giving 0
    return frac * float(np.sum(np.abs(inst.beta_true)))          # a fraction of ||beta*||_1


@pytest.mark.parametrize("kind,storage,restart", [(0, "f64", True), (1, "f64", True), (0, "f32", False),
                                                  (1, "f32", True)])
def test_lasso_trace_matches_oracle(dev, kind, storage, restart):
    import paper_2603_01306_amd as pr
    inst = make_instance(n=400, p=300, corr=0.7, k_true=8, snr=5.0, loss=0, seed=60 + kind, storage=storage)
    ctx = _ctx(dev, inst)
    lam = _lam(inst, kind, 0.1 if kind == 0 else 0.8)
    L = 2.02 * float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    its = 400
    tr = _trace(dev, its)
    method = pr.FISTA_GAP if restart else pr.FISTA
    r = ctx.lasso_solve(kind, lam, want_zeta=True, rel_gap_tol=1e-10, max_iter=its, L=L, method=method, trace=tr)
    ref = oracle.lasso_solve(inst.Xcm, inst.y, kind, lam, L=L, tol=1e-10, max_iter=its,
                             method=oracle.FISTA_GAP if restart else oracle.FISTA, trace_cap=its + 1)
    print({k: v for k, v in r.items() if k not in ("beta", "zeta")}, ref["iters"], ref["restarts"], flush=True)
    assert r["iters"] == ref["iters"] and r["restarts"] == ref["restarts"] and r["status"] == ref["status"]
    t = tr.cpu().numpy().reshape(-1, 2)[: r["iters"] + 1]
    scale = abs(ref["ub"])
    np.testing.assert_allclose(t[:, 0], ref["phi_trace"], rtol=0, atol=1e-10 * scale)
    np.testing.assert_allclose(t[:, 1], ref["phi_trace"] - ref["trace"], rtol=0, atol=1e-10 * scale)
    psi, s = oracle.lasso_dual(inst.Xcm, inst.y, kind, lam, r["zeta"].cpu().numpy())
    assert abs(psi - r["lower_bound"]) <= 1e-12 * scale and s == pytest.approx(1.0, abs=1e-12)
    b = r["beta"].cpu().numpy()
    phi = float(np.sum((inst.y - oracle.matvec(inst.Xcm, b)) ** 2)) + oracle.lasso_G(kind, b, lam)
    assert abs(phi - r["primal"]) <= 1e-12 * scale
    ctx.close()


@pytest.mark.parametrize("kind", [0, 1])
def test_lasso_full_size_certificate(dev, kind):
    """l1-regularised and l1-ball LASSO on the n = 16384, p = 8192 FP32 design
    to a 1e-6 gap with the gap restart: the oracle recomputes Psi at the
    returned dual point and Phi at the returned beta over the stored X."""
    import paper_2603_01306_amd as pr
    inst = config_instance("ls_root_n16384_p8192_f32")
    ctx = _ctx(dev, inst)
    lam = _lam(inst, kind, 0.05 if kind == 0 else 1.0)
    r = ctx.lasso_solve(kind, lam, want_zeta=True, max_iter=20000)
    print(kind, lam, {k: v for k, v in r.items() if k not in ("beta", "zeta")}, flush=True)
    assert r["status"] == pr.CONVERGED
    psi, _ = oracle.lasso_dual(inst.Xcm, inst.y, kind, lam, r["zeta"].cpu().numpy())
    b = r["beta"].cpu().numpy()
    phi = float(np.sum((inst.y - oracle.matvec(inst.Xcm, b)) ** 2)) + oracle.lasso_G(kind, b, lam)
    assert abs(psi - r["lower_bound"]) <= 1e-10 * abs(psi)
    assert abs(phi - r["primal"]) <= 1e-10 * abs(phi)
    assert 0.0 <= (phi - psi) / abs(phi) <= 1e-6
    ctx.close()


def test_lasso_rejects_bad_arguments(dev):
    import paper_2603_01306_amd as pr
    inst = make_instance(n=64, p=32, corr=0.5, k_true=3, snr=5.0, loss=1, seed=2, storage="f64")
    c = _ctx(dev, inst)
    with pytest.raises(pr.PrError):
        c.lasso_solve(pr.L1_REG, 1.0)                      # logistic context
    c.close()
    inst = make_instance(n=64, p=32, corr=0.5, k_true=3, snr=5.0, loss=0, seed=2, storage="f64")
    c = _ctx(dev, inst)
    for kind, lam, kw in ((2, 1.0, {}), (0, 0.0, {}), (0, 1.0, dict(method=pr.PGD))):
        with pytest.raises(pr.PrError):
            c.lasso_solve(kind, lam, **kw)
    c.close()
